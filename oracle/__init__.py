"""The oracle: a plain FP64 CPU reference tracker written from the paper.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import, load or run anything here.  It
shares no code with the GPU library.
"""
