"""MI355X-native occupancy-grid ray sampler: dense grid -> VDB tree ->
hierarchical DDA -> packed fixed-step samples, plus a fused volume-rendering
composite and a batched multi-scene launch.

Submodules: ``api`` (the Python binding of the C-ABI library, loaded on first
use) and ``scenes`` (seeded synthetic inputs).  Importing the package itself
touches no GPU and loads no library.
"""
