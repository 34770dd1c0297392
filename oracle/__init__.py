"""FP64 CPU oracle for the slice-streaming LJ path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``.  The product path never imports it.
"""
