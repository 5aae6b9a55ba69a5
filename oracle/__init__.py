"""Plain FP64 CPU oracle for the ADI-Newton thin-film step (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the GPU library.
"""
