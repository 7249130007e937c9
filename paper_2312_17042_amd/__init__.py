"""MI355X (gfx950) CTENO/CTENOZ finite-volume hot path: HIP kernels behind a C ABI.

Modules: ``cteno`` (ctypes binding of libcteno.so), ``workloads`` (seeded
synthetic meshes and exact solutions), ``build`` (hipcc build of the library).
"""
