"""SMMO (Single-Method Multiple-Objects) execution on AMD Instinct MI355X.

libsmmo.so (HIP, gfx950) implements the heap, the device allocator and the
do-all methods behind the C ABI in include/smmo.h; ``smmo`` is its Python
binding and ``sims`` drives the Game-of-Life, n-body and spring-mesh
workloads through it.
"""
