"""MI355X-native linear lattice Boltzmann acoustics (arXiv:1704.03172).

The compute path is the HIP library built from csrc/ (C-ABI declared in
include/lbwave.h); `lbwave` is its thin ctypes binding, with torch used only
for device memory and streams.  `inputs` builds seeded synthetic workloads.
Nothing is imported eagerly so that `inputs` can be used without a GPU.
"""
