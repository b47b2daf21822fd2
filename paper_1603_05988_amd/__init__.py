"""MI355X-native deflated Hutchinson / hierarchical-probing estimation of Tr(D^-1).

The computation lives in the HIP library libdhtrace.so (C ABI, include/dhtrace.h);
`paper_1603_05988_amd._lib` is its ctypes binding.  `workloads` generates the
seeded synthetic inputs.  Nothing here falls back to a CPU path: without the
built library the binding raises.
"""
__all__ = ["workloads"]
