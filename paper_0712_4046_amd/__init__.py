"""MI355X-native multipoint Kronecker substitution (exact products in Z[x] and (Z/pZ)[x]).

The product path is the HIP library libksmul.so (C ABI in include/ks.h); ``ks`` is its thin
Python binding and ``workloads`` draws seeded synthetic inputs.
"""
