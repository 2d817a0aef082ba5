"""SGF (sparse geometric factorization) preconditioned CG on AMD MI355X.

The compute path is the HIP library ``libsgf.so`` (C ABI in include/sgf.h);
``paper_1907_03406_amd.sgf`` is its ctypes binding.
"""
