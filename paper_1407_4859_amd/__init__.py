"""MI355X-native data-layout engine: layout remaps, layout-generic section
kernels and the two-level (per-section greedy, whole-program shortest path)
layout selection, behind the C-ABI library ``libadha.so``."""
