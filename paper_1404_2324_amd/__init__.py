"""MI355X-native hybrid symplectic N-body step (Grimm & Stadel, GENGA,
arXiv:1404.2324): hand-written gfx950 HIP kernels behind a C ABI
(``include/genga.h``), with a thin ctypes binding in ``genga``."""
