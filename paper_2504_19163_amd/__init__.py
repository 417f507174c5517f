"""Bernstein-bound caustics on AMD Instinct MI355X.

The method runs in the HIP library libbbc.so (C ABI in include/bbc.h); this
package holds its Python binding (bbc), its build step (build_lib) and the
seeded input generators (scenes).
"""
