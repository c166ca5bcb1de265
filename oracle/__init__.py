"""CPU oracle for batched Monte Carlo graph propagation (FS_GPlib, arxiv 2603.14895).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.

Two independent implementations of the same contract live here:

* ``fsg_oracle.c`` -- the plain loop nest of Algorithm 1 (per replicate, per
  step, per node, per in-edge) over uint8 states, plus a live-edge BFS for
  independent cascade; OpenMP over replicates only.  Wrapped by
  :mod:`oracle.native`.
* :mod:`oracle.twin` -- a pure-Python twin for tiny inputs (Philox on Python
  integers, dictionary-free list loops), used to cross-check the C code.

Pins that tie both to the paper and to mathematics (closed forms, exhaustive
enumeration of live-edge worlds, exact Markov chains, published Philox test
vectors) are in ``tests/test_oracle_*.py``.
"""
from . import native, twin  # noqa: F401
from .native import (  # noqa: F401
    IC, SI, SIS, SIR, LT, SEIR, SEIS, SWIR,
    IC_UNIFORM, IC_WEIGHTED_CASCADE, IC_PER_EDGE,
    DOM_IC_EDGE, DOM_NODE_STEP, DOM_LT_THRESH,
    philox4x32_10, draw, draw_many, thr, sir_table, simulate, ic_live_edge, hk, whk, hk_rows, build,
)
