"""MI355X-native batched acceptance-walk nested sampler (arXiv:2509.04336).

The compute path is the HIP library ``libnsmi.so`` behind the C ABI declared
in ``include/nsmi.h``; ``paper_2509_04336_amd.nsmi`` is its ctypes binding.
``paper_2509_04336_amd.inputs`` builds seeded synthetic workloads.
"""
__all__ = ["inputs", "nsmi"]
