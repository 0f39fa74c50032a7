"""MI355X-native FSMP: batched reversible-jump MCMC over PMT photo-electron sequences.

The sampler runs in hand-written HIP kernels for gfx950 behind the C ABI declared
in ``include/fsmp.h`` (``libfsmp.so``); :mod:`.fsmp` is a thin ctypes binding with
the same names.  :mod:`.synth` generates seeded synthetic workloads.
"""
