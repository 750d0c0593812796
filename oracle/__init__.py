"""CPU oracle for the ClusterMerge hot path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct implementations of
what the GPU library computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with ``paper_1908_10574_amd`` and never imports it.

Contents:
  * ``sw`` / ``sw_span`` / ``sw_batch`` / ``span_batch`` / ``traceback_batch``
    -- scalar Gotoh Smith-Waterman (score, end, start, alignment columns) in C
    (``sw_oracle.c``), loaded with ctypes;
  * ``brute`` -- enumeration of every local alignment (tiny inputs) and the
    cubic general-gap recurrence; used to pin the C code;
  * ``clustermerge`` -- Algorithm 1 (Cluster Set Merge) and Algorithm 2
    (BottomUpMerge) written out sequentially, the final in-cluster
    all-to-all and recall;
  * ``screen`` -- the hashed 3-mer featurizer and the MLP screen in numpy.
"""
from .sw import sw, sw_span, sw_batch, span_batch, traceback_batch, lib_path  # noqa: F401
