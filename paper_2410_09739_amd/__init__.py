"""MI355X-native D3Q27 Fokker-Planck central-moment lattice Boltzmann method.

The product is the C-ABI library ``liblbm.so`` (``include/lbm.h``), built from
``csrc/`` for gfx950.  ``paper_2410_09739_amd.lbm`` is its thin ctypes binding;
``paper_2410_09739_amd.workloads`` builds seeded synthetic inputs.  Submodules
are imported lazily so that importing the package touches no GPU.
"""
__all__ = ["lbm", "workloads"]
