"""CPU FP64 oracle for the periodic voxel homogenization path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it and shares no code with it; both sides only share the seeded
input generators of ``gmt_inputs``.

Everything here is plain numpy/scipy in float64, written from the paper's
definitions (Sec. 3.1 problem statement, Sec. 4.1 sparse hierarchy, Sec. 4.6
EBE operator and Galerkin coarse operators, Alg. 1/2 V-cycle, App. E transfer
operators, App. F homogenization).  Each module says which passage it follows.

Conventions fixed where the paper is silent:
* voxel arrays are indexed ``[z, y, x]``; linear index ``x + N*(y + N*z)``;
* active elements / nodes of a level are sorted by linear index, id = rank;
* hex8 local corner ``a + 2b + 4c`` sits at offset ``(a, b, c)``;
* DOF ``d`` of node ``i`` for load case ``m`` lives at ``u[i, m, d]``;
* Voigt order (11, 22, 33, 23, 13, 12) with engineering shear strains.

Parity status of each function is stated in its docstring; the network
reference (learned path) is the only part whose *quality* is parity unpinned.
"""
