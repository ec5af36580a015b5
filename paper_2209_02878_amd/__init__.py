"""MI355X-native (gfx950, HIP) segment / triangle-mesh intersection.

Tests N_r line segments against a triangle mesh through a linear BVH built on
the GPU, in three modes: a boolean crossing flag per segment, the first hit
(t, barycentric u and v, hit point, triangle id) and every crossing in a
bounded per-segment buffer with overflow retry.  The work runs in hand-written
HIP kernels behind a C ABI (include/rsi.h); `rsi` is the thin ctypes binding.
"""
