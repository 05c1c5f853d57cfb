"""MI355X-native Spring-Ising hot path (arXiv 2305.07187).

The compute lives in libspring_ising.so (hand-written HIP for gfx950) behind
the C ABI of include/spring_ising.h; ``spring_ising`` is its Python binding
and ``instances`` the seeded synthetic input generator.  Importing the
package does not load the library; the binding loads it on first use.
"""
__all__ = ["spring_ising", "instances", "build"]
