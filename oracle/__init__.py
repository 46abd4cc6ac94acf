"""The oracle: plain CPU references of what the GPU sorter computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import anything here; the product
path (``paper_1612_02557_amd``) never does, and shares no code with it.

* ``oracle_sort.c`` (C, built into ``liboracle.so``): stable LSD byte-wise
  counting sort (paper, Sec. 1), its T-thread form, one-digit histogram and
  one-digit stable partition, and duplicate removal with run counts over
  key-ordered records (the k-mer counting application, Sec. 5).
* ``mlp_ref`` (numpy, float64): the scheduler network's forward pass, loss,
  gradients and Adam step.
* ``sched_ref`` (Python): the heuristic procedure rules restated from the
  paper's thresholds (Sec. 3.2-3.5), and the regret of a choice.
* ``search_ref`` (Python): the suffix array of a text and the suffix-array
  range of each k-character query prefix (pattern search, Sec. 5).
"""
from .sort_ref import (  # noqa: F401
    lib,
    sort,
    sort_threads,
    sort_segments,
    partition,
    digit_histogram,
    count_runs,
    sort_count,
)
