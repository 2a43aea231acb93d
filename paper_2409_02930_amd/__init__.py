"""MI355X-native mean-field lattice Boltzmann for reactive mixtures in porous media.

The compute path is the HIP library built from ``csrc/`` (see ``build.py``);
``lbm`` is its ctypes binding.
"""
__all__ = ["lbm", "build"]
