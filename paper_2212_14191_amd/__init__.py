"""MI355X-native (gfx950) NTT / HMULT hot path of TensorFHE (arXiv 2212.14191).

The compute path is the C-ABI library ``libtfhe.so`` (hand-written HIP
kernels); ``paper_2212_14191_amd.tfhe`` is its thin ctypes binding.  Importing
the package itself loads nothing, so ``paper_2212_14191_amd.inputs`` (seeded
synthetic inputs) can be used without a GPU.
"""
