"""MI355X-native slice-streaming Lennard-Jones MD (cyclic data streaming, one GPU).

Importing the package loads nothing native; ``paper_2507_11289_amd.md`` binds the
HIP library and fails loudly when it is not built.
"""
__all__ = ["inputs"]
