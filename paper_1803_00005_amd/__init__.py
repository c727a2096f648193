"""MI355X-native hardware-efficient guided filter (HGF) for multi-label cost volumes.

``synth`` draws seeded synthetic workloads; ``hgf`` binds the HIP library
(``libhgf.so``, built by ``build_lib``) through its C ABI.
"""
__all__ = ["synth", "hgf", "build_lib"]
