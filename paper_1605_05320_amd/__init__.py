"""MI355X-native hot path of adjoint-guided refinement flagging for shallow-water
tsunami modelling: HIP kernels for gfx950 behind a C ABI (``include/swe.h``),
with a thin ctypes binding (``paper_1605_05320_amd.swe``)."""
