"""CPU FP64 oracle of the SGF factorization and SGF-preconditioned CG.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.
"""
