"""MI355X-native Blacklight hot path: camera, DP RK5(4) Kerr geodesics and
polarized thermal-synchrotron transfer in hand-written HIP kernels behind a
C ABI (libblgpu.so).  `blgpu` is the ctypes binding, `synth` the seeded input
generator."""
