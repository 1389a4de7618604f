"""CPU FP64 oracle for the PySchedCL attention / fork-join DAG path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this package: it is used by the
tests under ``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py``.  It shares no code with the HIP library (``paper_2009_07482_amd``); the two meet
only in the seeded input generators of ``workloads``, which hold none of the method's arithmetic.

Modules
  kernels    -- the four data-parallel kernels of the DAG in float64 (GEMM, transpose,
                row softmax, add), each the plain definition.
  bf16       -- round-to-nearest-even to bfloat16 and to float32, written from the IEEE /
                bfloat16 bit layouts.
  dag        -- executes a DAG spec in a topological order (Def. 5 of Sec. III); exact FP64 mode
                and a storage-dtype-emulating mode.
  attention  -- the multi-head attention layer of Sec. V written directly as formulas.
  validator  -- happens-before checker for exported command-queue structures (Def. 4, rules
                (i)-(iii) of Sec. III, Def. 5) and a brute-force interleaving checker.
  mlp        -- FP64 reference of the 3-layer MLP cost model: forward, MSE loss, backward,
                Adam.

Parity status: every function here is pinned by ``tests/test_oracle_*.py`` except the cost
model's makespan *predictions*, which have no published values (parity unpinned; they are assessed
by measured makespans instead).
"""
from . import kernels, bf16, dag, attention, validator, mlp  # noqa: F401
