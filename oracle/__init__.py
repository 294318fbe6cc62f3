"""Plain, slow FP64 CPU oracle of the two-level GenEO-type Schwarz method.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path may import, call or
link this package: only tests/, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP library; the only
common module is `workloads`, which generates the seeded inputs.

Every function cites the passage of Bootland, Dolean, Nataf & Tournier,
"A robust and adaptive GenEO-type domain decomposition preconditioner for
H(curl) problems in three-dimensional general topologies" (arXiv 2311.18783)
that it follows.  Where the method's result has a plain definition the
oracle writes that definition out with numpy / scipy primitives (dense
Cholesky, dense symmetric eigensolver, sparse LU); there is no blocking,
fusion or reordering beyond the definitions.

Pins (tests/test_oracle_*.py): K G = 0, element identities for constant and
linear fields, first-order convergence to a manufactured solution, the
paper's dof / NK / SNK counts (the SNK count through the overlapping
subdomains of Decomposition), hand-computed recursive-bisection parts,
overlap layers and smooth partition-of-unity values, the partition-of-unity
identity, k0 / k1 on geometries where they follow by hand, projector
identities, the GEVP bound lemma, the condition-number theorem (spectrum of
M^-1 A in [1/81, 8] on the 8^3 cube), brute-force dense cross-checks on tiny
meshes, GMRES against its defining minimal-residual property.  Parity
unpinned: none of the functions below; the MLP (oracle/mlp.py) has no
counterpart in the paper and is pinned by central finite differences.
"""
