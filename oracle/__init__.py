"""CPU oracle for the filtered Lanczos procedure: TEST INFRASTRUCTURE.

A plain FP64 implementation written from the paper.  Only ``tests/``, the
smoke check and the benchmark's CPU-baseline leg may use it; the GPU library
never imports, links or calls anything here.
"""
