"""MI355X-native matrix-free spectral-element PCG (FP64, mixed FP32/FP64,
iterative refinement, batched solves, learned flexible-CG preconditioner).

The compute path is the HIP library ``libmxsem.so`` behind the C ABI in
``include/mxsem.h``; ``paper_2503_02134_amd.mxsem`` is its Python binding.
Importing this package does not load the library; ``workloads`` (synthetic
inputs) is usable without a GPU.
"""
