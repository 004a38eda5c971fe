"""CPU oracle for the coupled point + field region grower.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(the HIP path) never imports, links or calls anything here, and nothing here
imports the product library: the two share only the seeded input generator.

Contents
  bfs    -- single-thread breadth-first grower in plain C (grow_bfs.c),
            loaded with ctypes; built by build_oracle().
  sweep  -- the fixed-point definition iterated literally: synchronous full
            sweeps F(X) = S_adm ∪ (Adm ∩ N(X)) in numpy until nothing changes.
  check  -- the invariants that single out the result, and an explicit edge
            list of the coupled graph for library connected-components.
  slic   -- the 4D clustering, cluster merging and feature statistics.
  segments -- the trajectory segment rule: runs of >= 2 consecutive steps
            of a particle in one feature.
"""
from .bfs import build_oracle, oracle_grow, oracle_grow_queries, oracle_seed_ids  # noqa: F401
from .sweep import sweep_grow  # noqa: F401
from .check import check_invariants, edge_list, components_grow, reach_grow  # noqa: F401
