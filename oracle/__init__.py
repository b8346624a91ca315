"""FP64 CPU oracle of the multilevel lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library
(no kernels, headers, tables or helpers); only the seeded input generators
in ``workloads`` feed both sides.

It is written to be plain and slow and to follow the paper step by step
(Qi, Klimach, Roller: "Implementation of the compact interpolation within
the octree based Lattice Boltzmann solver Musubi"):

* lattice.py  -- DdQq velocity sets and weights (Sec. 2.1)
* treeid.py   -- treeID decoding, Z-curve order, workload weights (Sec. 3.1)
* mesh.py     -- level-wise element lists, ghost classification, neighbour
                 and interpolation-source tables (Sec. 2.2, Sec. 3.2)
* physics.py  -- moments, equilibrium, strain rate, BGK (Sec. 2.1)
* interp.py   -- the four-source compact interpolation (Sec. 2.2,
                 Eqs. compact_3D_u / compact_3D_s, Steps 1-5)
* solver.py   -- recursive multilevel time stepping with NaN-poisoned
                 ghosts, diagnostics (Sec. 2.2, 2.3)
* tgv.py      -- Taylor-Green closed form and error norms (Sec. 4.1)
* adjoint.py  -- reverse pass of the whole oracle run by automatic
                 differentiation, plus central finite differences

Where the paper is silent or garbled, the reading taken is stated in the
docstring of the function that implements it.  Parity unpinned: the 2D
interpolation of non-quadratic data (the 2D algorithm is only referenced by
the paper), the choice of tetrahedron for non-quadratic data, the initial
ghost values and the far-field boundary conditions are fixed by those
readings alone.
"""
